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
//
// Direct mode (the default) copies nothing at stage time: the device keeps
// as many neighbour indices as the budget allows (a prefix of the CSR
// table), and the stage kernel reads the others across the host link from
// the pinned buffer itself, staging each workgroup's run of arcs in LDS with
// 16-byte loads.  One launch per stage, no copy stream, no events; measured
// on MI355X, such kernel reads of pinned memory move as many bytes per second
// as the copy engine (55 GB/s) and need no host work per tile.

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
  int mode = QW_STREAM_DIRECT;
  std::vector<int32_t> row;  // ring: tile t holds rows [row[t], row[t+1]); direct: workgroup tiles
  std::vector<int64_t> arc;  // ring: arcs [arc[t], arc[t+1])
  int64_t slot_arcs = 0;     // ring: neighbour indices per slot
  int64_t split = 0;         // direct: arcs [0, split) keep their indices on the device
  size_t rp_bytes = 0, bits_bytes = 0, mlist_bytes = 0, resident = 0, slot_stride = 0, wg_bytes = 0;
  size_t device_bytes = 0, host_bytes = 0;
};

int64_t round4(int64_t x) { return (x + 3) & ~int64_t{3}; }

// direct mode: workgroup tiles of at most kDirRows rows and kDirArcs arcs; a
// longer row is a tile of its own
void direct_tiles(const int32_t *rp, int64_t n, std::vector<int32_t> *row) {
  row->clear();
  int64_t r = 0;
  while (r < n) {
    row->push_back(static_cast<int32_t>(r));
    const int64_t r0 = r, a0 = rp[r];
    ++r;
    while (r < n && r - r0 < kDirRows && rp[r + 1] - a0 <= kDirArcs) ++r;
  }
  row->push_back(static_cast<int32_t>(n));
}

int schedule(const qw_plan *p, size_t budget, int mode, Schedule *out) {
  if (!p) return set_error(QW_EINVAL, "null plan");
  if (mode != QW_STREAM_DIRECT && mode != QW_STREAM_RING) return set_error(QW_EINVAL, "unknown stream mode %d", mode);
  if (p->kind != QW_CTQW || p->structure != kGeneral)
    return set_error(QW_EUNSUPPORTED, "out-of-core evolution needs a CTQW plan on the CSR path (QW_LAYOUT_CSR)");
  if (p->n == 0) return set_error(QW_EINVAL, "empty graph");
  Schedule &sc = *out;
  sc.mode = mode;
  sc.rp_bytes = sizeof(int32_t) * static_cast<size_t>(p->n + 1);
  sc.bits_bytes = sizeof(uint32_t) * static_cast<size_t>((p->n + 31) / 32);
  sc.mlist_bytes = sizeof(int32_t) * static_cast<size_t>(std::max<int32_t>(p->n_marked, 1));
  sc.resident = align256(sc.rp_bytes) + align256(sc.bits_bytes) + align256(sc.mlist_bytes);
  const size_t walk = p->state_bytes + p->work_bytes;
  const int32_t *rp = reinterpret_cast<const int32_t *>(p->image.data() + p->off_rp);
  if (mode == QW_STREAM_DIRECT) {
    direct_tiles(rp, p->n, &sc.row);
    sc.arc.clear();
    sc.wg_bytes = align256(sizeof(int32_t) * sc.row.size());
    const size_t fixed = walk + sc.resident + sc.wg_bytes;
    if (budget < fixed)
      return set_error(QW_ENOMEM,
                       "device budget of %zu bytes is below the state, workspace and resident tables (%zu bytes)",
                       budget, fixed);
    // the prefix takes whole 256-byte units of what is left (so the buffer stays
    // within the budget), or the whole padded table when that fits
    const int64_t padded = round4(p->n_arcs);
    const size_t left = budget - fixed;
    sc.split = align256(sizeof(int32_t) * static_cast<size_t>(padded)) <= left
                   ? padded
                   : static_cast<int64_t>((left & ~static_cast<size_t>(255)) / sizeof(int32_t));
    sc.device_bytes = sc.resident + sc.wg_bytes + align256(sizeof(int32_t) * static_cast<size_t>(sc.split));
    sc.host_bytes = sizeof(int32_t) * static_cast<size_t>(std::max<int64_t>(padded, 4));
    return QW_OK;
  }
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
  p->h_col_dev = nullptr;
  p->d_ring = nullptr;
  p->d_wg_row = nullptr;
  p->d_prefix = nullptr;
  p->st_n_wg = 0;
  p->st_split = 0;
}

int evolve_streamed(const qw_plan *p, void *psi, unsigned char *work, int64_t steps, double *d_p, double *d_norm,
                    double *d_pmarked, hipStream_t s) {
  const bool c128 = p->dtype == QW_C128;
  const GraphView &g = p->view;
  const int K = p->K;
  if (steps > 0 && p->st_mode == QW_STREAM_DIRECT) {
    void *w0 = work, *w1 = work + p->off_w1;
    for (int64_t i = 0; i < steps; ++i) {
      const void *yin = psi;
      for (int k = K; k >= 1; --k) {
        void *yout = (k == 1) ? (K == 1 ? w0 : psi) : (((K - k) & 1) ? w1 : w0);
        const double alpha = p->gamma * p->dt / k, beta = p->dt / k;
        QW_TRY(ctqw_direct_stage(c128, g, p->d_wg_row, p->st_n_wg, p->d_prefix, p->h_col_dev, p->st_split, yin, psi,
                                 yout, alpha, beta, s),
               "out-of-core CTQW stage kernel");
        yin = yout;
      }
      if (K == 1) QW_TRY(copy_state(c128, p->n, w0, psi, s), "state copy kernel");
    }
  } else if (steps > 0) {
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

int qw_plan_stream_sizes(const qw_plan *plan, size_t device_budget, int mode, size_t *host_bytes,
                         size_t *device_bytes, int64_t *n_tiles, int64_t *device_arcs) {
  Schedule sc;
  try {
    const int st = schedule(plan, device_budget, mode, &sc);
    if (st != QW_OK) return st;
  } catch (const std::bad_alloc &) {
    return set_error(QW_ENOMEM, "host allocation failed");
  }
  if (host_bytes) *host_bytes = sc.host_bytes;
  if (device_bytes) *device_bytes = sc.device_bytes;
  if (n_tiles) *n_tiles = static_cast<int64_t>(sc.row.size()) - 1;
  if (device_arcs) *device_arcs = mode == QW_STREAM_DIRECT ? std::min<int64_t>(sc.split, plan->n_arcs) : 0;
  return clear_error();
}

int qw_plan_upload_streamed(qw_plan *p, size_t device_budget, int mode, void *h_pinned, size_t host_bytes,
                            void *d_buf, size_t device_bytes, void *stream) {
  if (!p || !h_pinned || !d_buf) return set_error(QW_EINVAL, "null plan or buffer");
  Schedule sc;
  try {
    const int st = schedule(p, device_budget, mode, &sc);
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
  if (reinterpret_cast<uintptr_t>(h_pinned) % 16 != 0) return set_error(QW_EINVAL, "host buffer not 16-byte aligned");
  const int32_t *h_dev = nullptr;
  if (mode == QW_STREAM_DIRECT) {
    // the kernel reads the buffer itself: it must be pinned memory mapped for the device
    void *dp = nullptr;
    if (hipHostGetDevicePointer(&dp, h_pinned, 0) != hipSuccess || !dp) {
      (void)hipGetLastError();
      return set_error(QW_EINVAL, "host buffer is not pinned memory the device can read (hipHostMalloc)");
    }
    h_dev = static_cast<const int32_t *>(dp);
  }
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
  const size_t col_bytes = sizeof(int32_t) * static_cast<size_t>(p->n_arcs);
  std::memcpy(h_pinned, p->image.data() + p->off_col, col_bytes);
  std::memset(static_cast<unsigned char *>(h_pinned) + col_bytes, 0, sc.host_bytes - col_bytes);  // 16-byte tail
  if (mode == QW_STREAM_DIRECT) {
    const size_t o_wg = sc.resident, o_pre = sc.resident + sc.wg_bytes;
    QW_TRY(hipMemcpyAsync(base + o_wg, sc.row.data(), sizeof(int32_t) * sc.row.size(), hipMemcpyHostToDevice, s),
           "tile table upload");
    const size_t pre = sizeof(int32_t) * static_cast<size_t>(std::min<int64_t>(sc.split, p->n_arcs));
    if (pre > 0)
      QW_TRY(hipMemcpyAsync(base + o_pre, p->image.data() + p->off_col, pre, hipMemcpyHostToDevice, s),
             "neighbour prefix upload");
    if (sc.split > p->n_arcs)  // the prefix holds every arc: its 16-byte tail from the zeroed host tail
      QW_TRY(hipMemcpyAsync(base + o_pre + pre, static_cast<unsigned char *>(h_pinned) + col_bytes,
                            sizeof(int32_t) * static_cast<size_t>(sc.split) - pre, hipMemcpyHostToDevice, s),
             "neighbour prefix tail");
    p->d_wg_row = reinterpret_cast<int32_t *>(base + o_wg);
    p->st_n_wg = static_cast<int64_t>(sc.row.size()) - 1;
    p->d_prefix = reinterpret_cast<int32_t *>(base + o_pre);
    p->st_split = sc.split;
    p->h_col_dev = h_dev;
  } else {
    QW_TRY(hipStreamCreateWithFlags(&p->st_copy, hipStreamNonBlocking), "copy stream");
    p->st_free.assign(kSlots, nullptr);
    p->st_copied.assign(kSlots, nullptr);
    for (int i = 0; i < kSlots; ++i) {
      QW_TRY(hipEventCreateWithFlags(&p->st_free[i], hipEventDisableTiming), "ring event");
      QW_TRY(hipEventCreateWithFlags(&p->st_copied[i], hipEventDisableTiming), "ring event");
    }
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
  p->st_mode = mode;
  if (mode == QW_STREAM_RING) {
    p->st_row = std::move(sc.row);
    p->st_arc = std::move(sc.arc);
    p->st_slots = kSlots;
    p->st_slot_arcs = sc.slot_arcs;
    p->d_ring = reinterpret_cast<int32_t *>(base + sc.resident);
  } else {
    p->st_row.clear();
    p->st_arc.clear();
    p->st_slots = 0;
  }
  p->d_graph = base;
  p->streamed = true;
  return clear_error();
}

}  // extern "C"
