// qw_evolve_static: qw_evolve with the workspace taken from a device array of
// fixed size that this library holds, for callers that cannot allocate device
// memory.  The array is a file-scope __device__ symbol: each GPU the library
// runs on holds its own copy from module load until the process ends.  Host
// code never passes the symbol itself to a kernel (in host code its name is a
// host-side stand-in, not a device address); it asks the runtime for the
// address on each device once, with that device current, and passes that.

#include <mutex>

#include "qw_plan.h"
#include "qwalk.h"

namespace {

constexpr size_t kStaticScratchBytes = static_cast<size_t>(QW_STATIC_SCRATCH_BYTES);
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// This device's address of `scratch`, looked up on the device's first call.
int scratch_on(int dev, void **out) {
  if (dev < 0 || dev >= kMaxDevices) return qwk::set_error(QW_EDEVICE, "device %d out of range", dev);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    int cur = 0;
    hipError_t e = hipGetDevice(&cur);
    if (e == hipSuccess && cur != dev) e = hipSetDevice(dev);
    void *ptr = nullptr;
    if (e == hipSuccess) e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    const hipError_t back = (cur != dev) ? hipSetDevice(cur) : hipSuccess;
    if (e != hipSuccess)
      return qwk::set_error(QW_EDEVICE, "static scratch address on device %d: %s", dev, hipGetErrorString(e));
    if (back != hipSuccess)
      return qwk::set_error(QW_EDEVICE, "restoring device %d: %s", cur, hipGetErrorString(back));
    if (!ptr) return qwk::set_error(QW_EDEVICE, "static scratch on device %d has no address", dev);
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return QW_OK;
}

}  // namespace

extern "C" {

int qw_evolve_static(const qw_plan *p, void *d_psi, int64_t steps, double *d_p, double *d_norm, double *d_pmarked,
                     void *stream) {
  if (!p) return qwk::set_error(QW_EINVAL, "null plan");
  if (p->work_bytes > kStaticScratchBytes)
    return qwk::set_error(QW_ENOMEM,
                          "plan needs %zu bytes of workspace; the allocation-free entry point holds %zu "
                          "(QW_STATIC_SCRATCH_BYTES)",
                          p->work_bytes, kStaticScratchBytes);
  hipStream_t s = static_cast<hipStream_t>(stream);
  int dev = 0;
  const hipError_t e = s ? hipStreamGetDevice(s, &dev) : hipGetDevice(&dev);
  if (e != hipSuccess) return qwk::set_error(QW_EDEVICE, "device of the stream: %s", hipGetErrorString(e));
  void *work = nullptr;
  const int st = scratch_on(dev, &work);
  if (st != QW_OK) return st;
  return qw_evolve(p, d_psi, work, kStaticScratchBytes, steps, d_p, d_norm, d_pmarked, stream);
}

}  // extern "C"
