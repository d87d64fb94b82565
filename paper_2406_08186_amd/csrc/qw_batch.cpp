// Batched execution of many walks: the qw_batch_* half of the C ABI.
//
// A batch is a fixed table of slots.  Each launch of the batched kernel
// advances every active slot by one unit (a Horner stage of a CTQW step, or a
// coined step), so walks of very different sizes share launches and the
// per-launch work is the sum of theirs.  The launch sequence is captured once
// into a hipGraph and replayed; a device-side launch counter (advanced by the
// last workgroup of each launch) lets every replay find its place, and the
// host keeps a mirror of it.  Slots can be filled and emptied between runs
// (continuous batching); the host rebuilds the tile table, placing each
// walk's tiles on one XCD, and uploads the tables on the caller's stream.

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <numeric>
#include <vector>

#include "qw_internal.h"
#include "qw_plan.h"
#include "qwalk.h"

using namespace qwk;

namespace {

constexpr int kCoefStride = 128;  // doubles per slot: alpha[64], beta[64]
constexpr int kMaxGrid = 2048;    // 8 workgroups per CU at 256 CUs
constexpr int kLdsMaxGrid = 256;  // the LDS-staged kernel: one workgroup per CU (144-156 KiB of LDS each)
constexpr int kGraphChunk = 16;   // launches per captured graph

size_t align256(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }

struct ScheduleKey {
  int dtype;
  int64_t rows_bucket;
  int64_t deg_bucket;
  bool operator<(const ScheduleKey &o) const {
    return std::tie(dtype, rows_bucket, deg_bucket) < std::tie(o.dtype, o.rows_bucket, o.deg_bucket);
  }
};
struct Schedule {
  int rows, xcd, kernel;
};
std::mutex g_tune_mu;
std::map<ScheduleKey, Schedule> g_tune_cache;

}  // namespace

struct qw_batch {
  int32_t capacity = 0, max_tiles = 0, dtype = QW_C64;
  int32_t rows_per_tile = 1024;
  bool xcd_aware = true;
  int32_t stage_kernel = QW_BATCH_LDS;  // kernel for CTQW walks on the ELL layout of degree <= 8
  bool use_graph = true;  // qw_batch_run replays captured launches (else launches each directly)
  int grid = 8;      // workgroups of the gather kernel
  int grid_lds = 8;  // workgroups of the LDS-staged kernel
  // host staging
  std::vector<WalkSlot> slots;
  std::vector<const qw_plan *> plans;
  std::vector<int64_t> steps;
  std::vector<double> coefs;
  std::vector<TileEntry> table;   // tiles of the gather and structured kernels
  std::vector<TileEntry> ltable;  // tiles of the LDS-staged kernel
  int32_t n_tiles = 0, n_ltiles = 0;
  uint64_t L_host = 0;
  std::vector<char> needs_perm_in;  // structured coined slots staged since the last commit
  bool has_struct = false;          // any structured coined slot in the table (k_batch_struct runs)
  bool has_lds = false;             // any LDS-staged tile (k_batch_ell_lds runs, last in the unit)
  bool run_gather = true;           // k_batch_stage runs (it has tiles, or it advances the counter)
  // device binding
  unsigned char *d_buf = nullptr;
  size_t off_ctl = 0, off_slots = 0, off_coefs = 0, off_tiles = 0, off_ltiles = 0, off_ntiles = 0, bytes = 0;
  // pinned staging for table uploads, and the event that guards its reuse
  unsigned char *h_stage = nullptr;
  size_t stage_bytes = 0;
  hipEvent_t staged = nullptr;
  bool staged_pending = false;
  // graph replay
  hipStream_t capture = nullptr;
  hipGraphExec_t exec = nullptr;

  BatchCtl *ctl() const { return reinterpret_cast<BatchCtl *>(d_buf + off_ctl); }
  WalkSlot *dslots() const { return reinterpret_cast<WalkSlot *>(d_buf + off_slots); }
  double *dcoefs() const { return reinterpret_cast<double *>(d_buf + off_coefs); }
  TileEntry *dtiles() const { return reinterpret_cast<TileEntry *>(d_buf + off_tiles); }
  TileEntry *dltiles() const { return reinterpret_cast<TileEntry *>(d_buf + off_ltiles); }
  // tile counts: [0] the gather table, [1] the LDS-staged table
  int32_t *dntiles() const { return reinterpret_cast<int32_t *>(d_buf + off_ntiles); }
};

namespace {

int dev_fail(hipError_t e, const char *what) {
  return set_error(QW_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define QW_TRY(expr, what)                              \
  do {                                                  \
    hipError_t e_ = (expr);                             \
    if (e_ != hipSuccess) return dev_fail(e_, what);    \
  } while (0)

void layout(qw_batch *b) {
  size_t off = 0;
  auto sec = [&](size_t n) {
    const size_t o = off;
    off = align256(off + std::max<size_t>(n, 4));
    return o;
  };
  b->off_ctl = sec(sizeof(BatchCtl));
  b->off_slots = sec(sizeof(WalkSlot) * b->capacity);
  b->off_coefs = sec(sizeof(double) * kCoefStride * b->capacity);
  b->off_tiles = sec(sizeof(TileEntry) * b->max_tiles);
  b->off_ltiles = sec(sizeof(TileEntry) * b->max_tiles);
  b->off_ntiles = sec(2 * sizeof(int32_t));
  b->bytes = off;
}

// Host copy of a plan's coined tile boundaries (from its device image).
std::vector<int32_t> plan_tiles(const qw_plan *p) {
  std::vector<int32_t> t(static_cast<size_t>(p->n_tiles) + 1);
  std::memcpy(t.data(), p->image.data() + p->off_tiles, sizeof(int32_t) * t.size());
  return t;
}

std::vector<int32_t> plan_row_ptr(const qw_plan *p) {
  std::vector<int32_t> r(static_cast<size_t>(p->n) + 1);
  std::memcpy(r.data(), p->image.data() + p->off_rp, sizeof(int32_t) * r.size());
  return r;
}

int wait_stage(qw_batch *b) {
  if (b->staged_pending) {
    QW_TRY(hipEventSynchronize(b->staged), "batch staging wait");
    b->staged_pending = false;
  }
  return QW_OK;
}

// True when a slot's CTQW walk runs on the LDS-staged kernel.
bool lds_slot(const qw_batch *b, const WalkSlot &w) {
  // the LDS-staged kernel addresses the vector by 32-bit byte offsets and
  // stages it with 16-byte loads (aligned buffers, at least 16 bytes of state)
  const int64_t elem = b->dtype == QW_C128 ? 16 : 8;
  const bool aligned = ((reinterpret_cast<uintptr_t>(w.psi) | reinterpret_cast<uintptr_t>(w.w0) |
                         reinterpret_cast<uintptr_t>(w.w1)) & 15) == 0;
  return b->stage_kernel == QW_BATCH_LDS && w.kind == QW_CTQW && w.ell_d >= 1 && w.ell_d <= 8 &&
         static_cast<int64_t>(w.n) * elem < (int64_t{1} << 31) && static_cast<int64_t>(w.n) * elem >= 16 &&
         aligned;
}

// Lay out walks' tiles by XCD: longest walks first, each onto the XCD with
// the least load so far; entry 8 i + x is the i-th tile of XCD x's list, so a
// kernel whose grid is a multiple of 8 runs all of a walk's tiles on one XCD.
struct Item {
  int32_t slot;
  int64_t load;
  std::vector<TileEntry> tiles;
};
std::vector<TileEntry> lay_out(std::vector<Item> &items, bool xcd_aware) {
  std::vector<TileEntry> table;
  if (xcd_aware) {
    std::sort(items.begin(), items.end(), [](const Item &x, const Item &y) { return x.load > y.load; });
    std::vector<std::vector<TileEntry>> lists(8);
    int64_t load[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (const Item &it : items) {
      const int x = static_cast<int>(std::min_element(load, load + 8) - load);
      load[x] += it.load;
      lists[x].insert(lists[x].end(), it.tiles.begin(), it.tiles.end());
    }
    size_t m = 0;
    for (const auto &l : lists) m = std::max(m, l.size());
    table.assign(8 * m, TileEntry{-1, 0, 0, 0});
    for (int x = 0; x < 8; ++x)
      for (size_t i = 0; i < lists[x].size(); ++i) table[8 * i + x] = lists[x][i];
  } else {
    for (const Item &it : items) table.insert(table.end(), it.tiles.begin(), it.tiles.end());
  }
  return table;
}

// Rebuild the tile tables from the active slots.
int build_table(qw_batch *b) {
  std::vector<Item> items, litems;
  for (int s = 0; s < b->capacity; ++s) {
    const WalkSlot &w = b->slots[s];
    if (w.kind < 0) continue;
    Item it;
    it.slot = s;
    const qw_plan *p = b->plans[s];
    if (w.kind == QW_CTQW) {
      const bool lds = lds_slot(b, w);
      const int R = lds ? (b->dtype == QW_C128 ? kLdsTileRows128 : kLdsTileRows64) : b->rows_per_tile;
      for (int64_t r = 0; r < p->n; r += R)
        it.tiles.push_back({s, static_cast<int32_t>(r), static_cast<int32_t>(std::min<int64_t>(p->n, r + R)), 0});
      it.load = p->n_arcs + 3 * p->n;
      if (lds) {
        litems.push_back(std::move(it));
        continue;
      }
    } else if (w.structure != kGeneral) {
      const int R = b->rows_per_tile;
      for (int64_t v = 0; v < p->n; v += R)
        it.tiles.push_back({s, static_cast<int32_t>(v), static_cast<int32_t>(std::min<int64_t>(p->n, v + R)), 0});
      it.load = 2 * p->n_arcs;
    } else {
      const std::vector<int32_t> t = plan_tiles(p);
      for (int32_t i = 0; i + 1 < static_cast<int32_t>(t.size()); ++i) it.tiles.push_back({s, t[i], t[i + 1], 0});
      it.load = 2 * p->n_arcs;
    }
    items.push_back(std::move(it));
  }
  bool has_struct = false;
  for (int s = 0; s < b->capacity; ++s)
    has_struct |= b->slots[s].kind == QW_COINED && b->slots[s].structure != kGeneral;
  std::vector<TileEntry> table = lay_out(items, b->xcd_aware);
  std::vector<TileEntry> ltable = lay_out(litems, b->xcd_aware);
  if (static_cast<int64_t>(table.size()) > b->max_tiles || static_cast<int64_t>(ltable.size()) > b->max_tiles)
    return set_error(QW_ENOMEM, "batch needs %zu + %zu tiles, capacity is %d per table", table.size(),
                     ltable.size(), b->max_tiles);
  const bool has_lds = !ltable.empty();
  // k_batch_stage runs when it has tiles, and also when nothing else would
  // advance the launch counter
  const bool run_gather = !table.empty() || !has_lds;
  // grids: multiples of 8 (keeps the XCD placement), no larger than the work
  const int grid = std::max(8, std::min(kMaxGrid, (static_cast<int>(table.size()) + 7) / 8 * 8));
  const int grid_lds = std::max(8, std::min(kLdsMaxGrid, (static_cast<int>(ltable.size()) + 7) / 8 * 8));
  if (has_struct != b->has_struct || has_lds != b->has_lds || run_gather != b->run_gather || grid != b->grid ||
      grid_lds != b->grid_lds) {
    if (b->exec) {
      (void)hipGraphExecDestroy(b->exec);  // the launch unit changed: re-captured at the next run
      b->exec = nullptr;
    }
  }
  b->has_struct = has_struct;
  b->has_lds = has_lds;
  b->run_gather = run_gather;
  b->grid = grid;
  b->grid_lds = grid_lds;
  b->table = std::move(table);
  b->ltable = std::move(ltable);
  b->n_tiles = static_cast<int32_t>(b->table.size());
  b->n_ltiles = static_cast<int32_t>(b->ltable.size());
  return QW_OK;
}

int upload_tables(qw_batch *b, hipStream_t s) {
  int st = wait_stage(b);
  if (st != QW_OK) return st;
  const size_t sl = sizeof(WalkSlot) * b->capacity;
  const size_t co = sizeof(double) * kCoefStride * b->capacity;
  const size_t ti = sizeof(TileEntry) * b->table.size();
  const size_t lt = sizeof(TileEntry) * b->ltable.size();
  unsigned char *h = b->h_stage;
  const size_t o_cnt = sl + co, o_ti = o_cnt + 256, o_lt = align256(o_ti + ti);
  std::memcpy(h, b->slots.data(), sl);
  std::memcpy(h + sl, b->coefs.data(), co);
  const int32_t counts[2] = {b->n_tiles, b->n_ltiles};
  std::memcpy(h + o_cnt, counts, sizeof counts);
  if (ti) std::memcpy(h + o_ti, b->table.data(), ti);
  if (lt) std::memcpy(h + o_lt, b->ltable.data(), lt);
  QW_TRY(hipMemcpyAsync(b->dslots(), h, sl, hipMemcpyHostToDevice, s), "batch slot upload");
  QW_TRY(hipMemcpyAsync(b->dcoefs(), h + sl, co, hipMemcpyHostToDevice, s), "batch coefficient upload");
  QW_TRY(hipMemcpyAsync(b->dntiles(), h + o_cnt, sizeof counts, hipMemcpyHostToDevice, s), "batch count upload");
  if (ti) QW_TRY(hipMemcpyAsync(b->dtiles(), h + o_ti, ti, hipMemcpyHostToDevice, s), "batch tile upload");
  if (lt) QW_TRY(hipMemcpyAsync(b->dltiles(), h + o_lt, lt, hipMemcpyHostToDevice, s), "batch tile upload");
  QW_TRY(hipEventRecord(b->staged, s), "batch staging event");
  b->staged_pending = true;
  return QW_OK;
}

int set_probe(qw_batch *b, unsigned int on, hipStream_t s) {
  int st = wait_stage(b);
  if (st != QW_OK) return st;
  std::memcpy(b->h_stage, &on, sizeof on);
  QW_TRY(hipMemcpyAsync(reinterpret_cast<unsigned char *>(b->ctl()) + offsetof(BatchCtl, probe), b->h_stage,
                        sizeof on, hipMemcpyHostToDevice, s),
         "batch probe flag");
  QW_TRY(hipEventRecord(b->staged, s), "batch staging event");
  b->staged_pending = true;
  return QW_OK;
}

// One batched unit: the structured coined tiles, then the gather kernel's
// tiles, then the LDS-staged tiles; the last kernel of the unit advances the
// launch counter.
hipError_t launch_one(qw_batch *b, hipStream_t s) {
  const bool c128 = b->dtype == QW_C128;
  if (b->has_struct) {
    const hipError_t e = batch_struct(c128, b->ctl(), b->dslots(), b->dtiles(), b->dntiles(), b->grid, s);
    if (e != hipSuccess) return e;
  }
  if (b->run_gather) {
    const hipError_t e =
        batch_stage(c128, b->ctl(), b->dslots(), b->dtiles(), b->dntiles(), b->grid, b->has_lds ? 0 : 1, s);
    if (e != hipSuccess) return e;
  }
  if (b->has_lds) return batch_ell_lds(c128, b->ctl(), b->dslots(), b->dltiles(), b->dntiles() + 1, b->grid_lds, 1, s);
  return hipSuccess;
}

int check_batch(const qw_batch *b) {
  if (!b) return set_error(QW_EINVAL, "null batch");
  if (!b->d_buf) return set_error(QW_ESTATE, "batch not bound (call qw_batch_bind first)");
  return QW_OK;
}

}  // namespace

extern "C" {

int qw_batch_create(int32_t capacity, int32_t max_tiles, int32_t dtype, qw_batch **out) {
  if (!out) return set_error(QW_EINVAL, "null output pointer");
  *out = nullptr;
  if (capacity < 1 || capacity > (1 << 20)) return set_error(QW_EINVAL, "capacity %d out of range", capacity);
  if (max_tiles < 8 || max_tiles > (1 << 28)) return set_error(QW_EINVAL, "max_tiles %d out of range", max_tiles);
  if (dtype != QW_C64 && dtype != QW_C128) return set_error(QW_EINVAL, "bad dtype %d", dtype);
  try {
    auto *b = new qw_batch();
    b->capacity = capacity;
    b->max_tiles = (max_tiles + 7) / 8 * 8;
    b->dtype = dtype;
    b->slots.assign(capacity, WalkSlot());
    for (auto &w : b->slots) w.kind = -1;
    b->plans.assign(capacity, nullptr);
    b->steps.assign(capacity, 0);
    b->needs_perm_in.assign(capacity, 0);
    b->coefs.assign(static_cast<size_t>(capacity) * kCoefStride, 0.0);
    b->grid = std::min(kMaxGrid, b->max_tiles);
    layout(b);
    *out = b;
  } catch (const std::bad_alloc &) {
    return set_error(QW_ENOMEM, "host allocation failed");
  }
  return clear_error();
}

int qw_batch_destroy(qw_batch *b) {
  if (!b) return clear_error();
  if (b->staged_pending) (void)hipEventSynchronize(b->staged);
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->capture) (void)hipStreamDestroy(b->capture);
  if (b->staged) (void)hipEventDestroy(b->staged);
  if (b->h_stage) (void)hipHostFree(b->h_stage);
  delete b;
  return clear_error();
}

int qw_batch_device_bytes(const qw_batch *b, size_t *bytes) {
  if (!b || !bytes) return set_error(QW_EINVAL, "null argument");
  *bytes = b->bytes;
  return clear_error();
}

int qw_batch_bind(qw_batch *b, void *d_buf, size_t bytes, void *stream) {
  if (!b || !d_buf) return set_error(QW_EINVAL, "null batch or buffer");
  if (bytes < b->bytes) return set_error(QW_ENOMEM, "batch buffer of %zu bytes, needs %zu", bytes, b->bytes);
  if (reinterpret_cast<uintptr_t>(d_buf) % 256) return set_error(QW_EINVAL, "batch buffer not 256-byte aligned");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (!b->h_stage) {
    b->stage_bytes = sizeof(WalkSlot) * b->capacity + sizeof(double) * kCoefStride * b->capacity + 256 +
                     2 * (sizeof(TileEntry) * b->max_tiles + 256) + 256;
    QW_TRY(hipHostMalloc(reinterpret_cast<void **>(&b->h_stage), b->stage_bytes, hipHostMallocDefault),
           "pinned staging allocation");
    QW_TRY(hipEventCreateWithFlags(&b->staged, hipEventDisableTiming), "batch event");
    QW_TRY(hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking), "batch capture stream");
  }
  if (b->exec) {
    (void)hipGraphExecDestroy(b->exec);
    b->exec = nullptr;
  }
  b->d_buf = static_cast<unsigned char *>(d_buf);
  int st = wait_stage(b);
  if (st != QW_OK) return st;
  BatchCtl zero{};
  std::memcpy(b->h_stage + b->stage_bytes - 256, &zero, sizeof zero);
  QW_TRY(hipMemcpyAsync(b->ctl(), b->h_stage + b->stage_bytes - 256, sizeof zero, hipMemcpyHostToDevice, s),
         "batch control reset");
  b->L_host = 0;
  for (int i = 0; i < b->capacity; ++i) {
    b->slots[i] = WalkSlot();
    b->slots[i].kind = -1;
    b->plans[i] = nullptr;
  }
  b->table.clear();
  b->ltable.clear();
  b->n_tiles = b->n_ltiles = 0;
  st = upload_tables(b, s);
  return st == QW_OK ? clear_error() : st;
}

int qw_batch_set_slot(qw_batch *b, int32_t slot, const qw_plan *p, void *d_psi, void *d_work,
                      size_t work_bytes, int64_t steps, double *d_hist) {
  int st = check_batch(b);
  if (st != QW_OK) return st;
  if (slot < 0 || slot >= b->capacity) return set_error(QW_EINVAL, "slot %d out of range", slot);
  if (!p || !d_psi || !d_work) return set_error(QW_EINVAL, "null plan, state or workspace");
  if (!p->d_graph) return set_error(QW_ESTATE, "plan not uploaded");
  if (p->streamed) return set_error(QW_EUNSUPPORTED, "plans bound for out-of-core evolution cannot join a batch");
  if (p->dtype != b->dtype) return set_error(QW_EINVAL, "plan dtype differs from the batch's");
  if (p->kind == QW_STAGGERED) return set_error(QW_EUNSUPPORTED, "staggered walks cannot join a batch");
  const bool coined_struct = p->kind == QW_COINED &&
                             (p->structure == kCycle || p->structure == kTorus || p->structure == kHypercube);
  if (!(p->structure == kGeneral || (p->kind == QW_CTQW && p->structure == kEll) || coined_struct))
    return set_error(QW_EUNSUPPORTED,
                     "batched walks need CSR plans, CTQW plans on the ELL path, or coined plans on a "
                     "cycle, torus or hypercube path");
  if (p->lattice() || p->coin == QW_SZEGEDY)
    return set_error(QW_EUNSUPPORTED,
                     "Fourier, matrix and Szegedy coins and the persistent shift cannot join a batch");
  if (work_bytes < p->work_bytes) return set_error(QW_ENOMEM, "workspace too small for the plan");
  if (steps < 0) return set_error(QW_EINVAL, "negative steps");
  if (p->n == 0) return set_error(QW_EINVAL, "empty graph");
  WalkSlot w;
  w.kind = p->kind;
  w.n = static_cast<int32_t>(p->n);
  w.K = p->kind == QW_CTQW ? p->K : 1;
  w.hadamard = p->coin == QW_HADAMARD;
  w.L0 = static_cast<int64_t>(b->L_host);
  w.units = steps * w.K;
  w.rp = p->view.rp;
  w.col = p->view.col;
  w.ell_d = p->structure == kEll ? p->view.ell_d : 0;
  w.pad0 = 0;
  w.structure = coined_struct ? p->structure : kGeneral;
  w.sdims[0] = p->dims[0];
  w.sdims[1] = p->dims[1];
  w.pad1 = 0;
  w.rev = p->view.rev;
  w.markbits = p->view.markbits;
  w.psi = d_psi;
  w.w0 = d_work;
  w.w1 = static_cast<unsigned char *>(d_work) + p->off_w1;
  w.hist = nullptr;
  double *co = b->coefs.data() + static_cast<size_t>(slot) * kCoefStride;
  std::fill(co, co + kCoefStride, 0.0);
  if (p->kind == QW_CTQW) {
    if (p->K < 2) return set_error(QW_EUNSUPPORTED, "batched CTQW needs Taylor order >= 2");
    for (int k = 1; k <= p->K; ++k) {
      co[k - 1] = p->gamma * p->dt / k;
      co[64 + k - 1] = p->dt / k;
    }
    w.hist = d_hist;
  } else {
    const std::vector<int32_t> t = plan_tiles(p);
    const std::vector<int32_t> rp = plan_row_ptr(p);
    for (size_t i = 0; i + 1 < t.size(); ++i)
      if (rp[t[i + 1]] - rp[t[i]] > kTileArcs)
        return set_error(QW_EUNSUPPORTED, "batched coined walks need every vertex degree <= %d", kTileArcs);
  }
  if (b->d_buf) {
    w.alpha = b->dcoefs() + static_cast<size_t>(slot) * kCoefStride;
    w.beta = w.alpha + 64;
  }
  b->slots[slot] = w;
  b->plans[slot] = p;
  b->steps[slot] = steps;
  b->needs_perm_in[slot] = coined_struct;
  return clear_error();
}

int qw_batch_clear_slot(qw_batch *b, int32_t slot) {
  if (!b) return set_error(QW_EINVAL, "null batch");
  if (slot < 0 || slot >= b->capacity) return set_error(QW_EINVAL, "slot %d out of range", slot);
  b->slots[slot] = WalkSlot();
  b->slots[slot].kind = -1;
  b->plans[slot] = nullptr;
  b->steps[slot] = 0;
  b->needs_perm_in[slot] = 0;
  return clear_error();
}

int qw_batch_commit(qw_batch *b, void *stream) {
  int st = check_batch(b);
  if (st != QW_OK) return st;
  st = build_table(b);
  if (st != QW_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  for (int i = 0; i < b->capacity; ++i) {
    if (!b->needs_perm_in[i]) continue;
    const qw_plan *p = b->plans[i];
    QW_TRY(coined_perm_in(b->dtype == QW_C128, p->view, b->slots[i].psi, b->slots[i].w0, s),
           "layout permutation kernel");
    b->needs_perm_in[i] = 0;
  }
  st = upload_tables(b, s);
  return st == QW_OK ? clear_error() : st;
}

int qw_batch_run(qw_batch *b, int64_t launches, void *stream) {
  int st = check_batch(b);
  if (st != QW_OK) return st;
  if (launches < 0) return set_error(QW_EINVAL, "negative launch count");
  hipStream_t s = static_cast<hipStream_t>(stream);
  int64_t replays = 0, direct = 0;
  qw_batch_launch_plan(b, launches, &replays, &direct);
  if (replays > 0) {
    if (!b->exec) {
      hipGraph_t g = nullptr;
      QW_TRY(hipStreamBeginCapture(b->capture, hipStreamCaptureModeRelaxed), "batch graph capture begin");
      hipError_t le = hipSuccess;
      for (int i = 0; i < kGraphChunk && le == hipSuccess; ++i) le = launch_one(b, b->capture);
      hipError_t ce = hipStreamEndCapture(b->capture, &g);
      if (le != hipSuccess) return dev_fail(le, "batch graph capture launch");
      if (ce != hipSuccess) return dev_fail(ce, "batch graph capture end");
      hipError_t ie = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (ie != hipSuccess) {
        b->exec = nullptr;
        return dev_fail(ie, "batch graph instantiate");
      }
    }
    for (int64_t i = 0; i < replays; ++i) QW_TRY(hipGraphLaunch(b->exec, s), "batch graph launch");
  }
  for (int64_t i = 0; i < direct; ++i) QW_TRY(launch_one(b, s), "batched stage kernel");
  b->L_host += static_cast<uint64_t>(launches);
  return clear_error();
}

int qw_batch_set_replay(qw_batch *b, int32_t use_graph) {
  if (!b) return set_error(QW_EINVAL, "null batch");
  b->use_graph = use_graph != 0;
  return clear_error();
}

int qw_batch_launch_plan(const qw_batch *b, int64_t launches, int64_t *graph_replays, int64_t *direct_launches) {
  if (!b) return set_error(QW_EINVAL, "null batch");
  if (launches < 0) return set_error(QW_EINVAL, "negative launch count");
  const int64_t replays = b->use_graph ? launches / kGraphChunk : 0;
  if (graph_replays) *graph_replays = replays;
  if (direct_launches) *direct_launches = launches - replays * kGraphChunk;
  return clear_error();
}

int qw_batch_remaining(const qw_batch *b, int32_t slot, int64_t *remaining) {
  if (!b || !remaining) return set_error(QW_EINVAL, "null argument");
  if (slot < 0 || slot >= b->capacity) return set_error(QW_EINVAL, "slot %d out of range", slot);
  const WalkSlot &w = b->slots[slot];
  if (w.kind < 0) {
    *remaining = 0;
  } else {
    const int64_t done = static_cast<int64_t>(b->L_host) - w.L0;
    *remaining = std::max<int64_t>(0, w.units - done);
  }
  return clear_error();
}

int qw_batch_launches(const qw_batch *b, int64_t *launches) {
  if (!b || !launches) return set_error(QW_EINVAL, "null argument");
  *launches = static_cast<int64_t>(b->L_host);
  return clear_error();
}

int qw_batch_readout(qw_batch *b, int32_t slot, double *d_p, double *d_norm, double *d_pmarked, void *stream) {
  int st = check_batch(b);
  if (st != QW_OK) return st;
  if (slot < 0 || slot >= b->capacity || b->slots[slot].kind < 0)
    return set_error(QW_EINVAL, "slot %d is empty or out of range", slot);
  int64_t rem = 0;
  qw_batch_remaining(b, slot, &rem);
  if (rem != 0) return set_error(QW_ESTATE, "slot %d still has %lld launches to run", slot, (long long)rem);
  const WalkSlot &w = b->slots[slot];
  const qw_plan *p = b->plans[slot];
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (w.kind == QW_COINED && w.structure != kGeneral) {
    // slot-major state: units alternate w0 -> w1 -> w0, so it ends in w1 after an odd count
    const void *fin = (b->steps[slot] & 1) ? w.w1 : w.w0;
    st = plan_struct_out(p, fin, w.psi, static_cast<unsigned char *>(w.w0), d_p, d_norm, d_pmarked, s);
    return st == QW_OK ? clear_error() : st;
  }
  if (w.kind == QW_COINED && (b->steps[slot] & 1))
    QW_TRY(copy_state(b->dtype == QW_C128, p->n_arcs, w.w0, w.psi, s), "state copy kernel");
  st = plan_readout(p, w.psi, static_cast<unsigned char *>(w.w0), d_p, d_norm, d_pmarked, s);
  return st == QW_OK ? clear_error() : st;
}

int qw_batch_set_schedule(qw_batch *b, int32_t rows_per_tile, int32_t xcd_aware) {
  if (!b) return set_error(QW_EINVAL, "null batch");
  if (rows_per_tile < 64 || rows_per_tile > (1 << 20)) return set_error(QW_EINVAL, "rows_per_tile out of range");
  b->rows_per_tile = rows_per_tile;
  b->xcd_aware = xcd_aware != 0;
  return clear_error();
}

int qw_batch_set_stage_kernel(qw_batch *b, int32_t kernel) {
  if (!b) return set_error(QW_EINVAL, "null batch");
  if (kernel != QW_BATCH_GATHER && kernel != QW_BATCH_LDS) return set_error(QW_EINVAL, "bad stage kernel %d", kernel);
  b->stage_kernel = kernel;
  return clear_error();
}

int qw_batch_get_schedule(const qw_batch *b, int32_t *rows_per_tile, int32_t *xcd_aware, int32_t *kernel) {
  if (!b) return set_error(QW_EINVAL, "null batch");
  if (rows_per_tile) *rows_per_tile = b->rows_per_tile;
  if (xcd_aware) *xcd_aware = b->xcd_aware;
  if (kernel) *kernel = b->stage_kernel;
  return clear_error();
}

int qw_batch_autotune(qw_batch *b, int32_t reps, void *stream, int32_t *rows_per_tile, int32_t *xcd_aware,
                      double *ms_per_launch) {
  int st = check_batch(b);
  if (st != QW_OK) return st;
  if (reps < 1) return set_error(QW_EINVAL, "reps must be >= 1");
  int64_t rows = 0, arcs = 0, walks = 0;
  bool any_ell8 = false, any_other = false;
  for (int s = 0; s < b->capacity; ++s) {
    const WalkSlot &w = b->slots[s];
    if (w.kind < 0) continue;
    if (b->L_host != static_cast<uint64_t>(w.L0))
      return set_error(QW_ESTATE, "autotune needs every active walk at its first unit (slot %d has started)", s);
    rows += b->plans[s]->n;
    arcs += b->plans[s]->n_arcs;
    ++walks;
    const bool ell8 = w.kind == QW_CTQW && w.ell_d >= 1 && w.ell_d <= 8;
    any_ell8 |= ell8;
    any_other |= !ell8;
  }
  if (walks == 0) return set_error(QW_ESTATE, "no active walks to tune on");
  const ScheduleKey key{b->dtype, static_cast<int64_t>(std::log2(static_cast<double>(rows))),
                        static_cast<int64_t>(std::lround(2.0 * arcs / rows))};
  hipStream_t s = static_cast<hipStream_t>(stream);
  auto finish = [&](double ms) {
    if (rows_per_tile) *rows_per_tile = b->rows_per_tile;
    if (xcd_aware) *xcd_aware = b->xcd_aware;
    if (ms_per_launch) *ms_per_launch = ms;
    int r = build_table(b);
    if (r == QW_OK) r = upload_tables(b, s);
    return r == QW_OK ? clear_error() : r;
  };
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end()) {
      b->rows_per_tile = it->second.rows;
      b->xcd_aware = it->second.xcd != 0;
      b->stage_kernel = it->second.kernel;
      return finish(-1.0);
    }
  }
  hipEvent_t e0, e1;
  QW_TRY(hipEventCreate(&e0), "event");
  QW_TRY(hipEventCreate(&e1), "event");
  st = set_probe(b, 1u, s);
  double best = 1e300;
  Schedule bestc{b->rows_per_tile, b->xcd_aware, b->stage_kernel};
  const int cand_r[] = {256, 512, 1024, 2048, 4096};
  const int cand_k[] = {QW_BATCH_LDS, QW_BATCH_GATHER};
  for (int kern : cand_k) {
    if (kern == QW_BATCH_LDS && !any_ell8) continue;  // the same schedules as the gather kernel
    for (int xi = 1; xi >= 0 && st == QW_OK; --xi) {
      for (int r : cand_r) {
        // with every walk on the LDS-staged kernel, rows per tile change nothing
        if (kern == QW_BATCH_LDS && !any_other && r != cand_r[0]) continue;
        b->rows_per_tile = r;
        b->xcd_aware = xi != 0;
        b->stage_kernel = kern;
        st = build_table(b);
        if (st == QW_ENOMEM) {  // this schedule's tile table does not fit max_tiles: skip it
          st = QW_OK;
          continue;
        }
        if (st == QW_OK) st = upload_tables(b, s);
        if (st != QW_OK) break;
        hipError_t e = launch_one(b, s);
        if (e == hipSuccess) e = hipEventRecord(e0, s);
        for (int i = 0; i < reps && e == hipSuccess; ++i) e = launch_one(b, s);
        if (e == hipSuccess) e = hipEventRecord(e1, s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) {
          st = dev_fail(e, "autotune probe");
          break;
        }
        const double per = ms / reps;
        if (per < best) {
          best = per;
          bestc = {r, xi, kern};
        }
      }
    }
  }
  const int st2 = set_probe(b, 0u, s);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != QW_OK) return st;
  if (st2 != QW_OK) return st2;
  if (best > 1e299) return set_error(QW_ENOMEM, "no candidate schedule fits max_tiles");
  b->rows_per_tile = bestc.rows;
  b->xcd_aware = bestc.xcd != 0;
  b->stage_kernel = bestc.kernel;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[key] = bestc;
  }
  return finish(best);
}

}  // extern "C"
