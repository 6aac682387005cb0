// noalloc.hip -- phgrms_denoise_noalloc: the pass loop of
// phgrms_denoise_async with its workspace in a fixed device array of the
// library, for callers that cannot allocate device memory (code under graph
// capture, tight serving loops, harnesses that forbid allocation).
//
// The array is a file-scope __device__ symbol: each GPU the library runs
// on holds its own copy until the process ends.  In host code its name is
// only a host-side stand-in, so the device address is looked up once per
// device with hipGetSymbolAddress and used everywhere instead.
#include <hip/hip_runtime.h>

#include <mutex>

#include "phgrms.h"
#include "phgrms_internal.hpp"

namespace {

static __device__ __align__(256) uint8_t scratch[PHGRMS_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on the current device (looked up on the
// first call there).
int scratch_address(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return phg::hip_fail(e, "current device");
  if (dev < 0 || dev >= kMaxDevices)
    return phg::fail(PHGRMS_EUNSUPPORTED, "device %d beyond the %d the library tracks", dev, kMaxDevices);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return phg::hip_fail(e, "scratch symbol address");
    if (p == nullptr) return phg::fail(PHGRMS_EDEVICE, "scratch symbol has no device address");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return PHGRMS_OK;
}

}  // namespace

extern "C" int phgrms_denoise_noalloc(const uint8_t* d_in, uint8_t* d_out, phgrms_params p,
                                      int64_t* d_changed, int32_t* d_iterations, void* stream) {
  int rc = phg::validate_params(p);
  if (rc != PHGRMS_OK) return rc;
  const phg::WsLayout l = phg::ws_layout(p);
  if (l.total > size_t(PHGRMS_NOALLOC_SCRATCH_BYTES))
    return phg::fail(PHGRMS_ENOSPC,
                     "a %dx%d image with k = %d needs %zu bytes of workspace; the library's fixed "
                     "scratch holds %zu (use phgrms_denoise_async with a workspace)",
                     p.rows, p.cols, p.k, l.total, size_t(PHGRMS_NOALLOC_SCRATCH_BYTES));
  void* ws = nullptr;
  if ((rc = scratch_address(&ws)) != PHGRMS_OK) return rc;
  // the same path as phgrms_denoise_async, over the fixed scratch (which
  // the pass loop clears where it must start at zero)
  return phgrms_denoise_async(d_in, d_out, p, ws, size_t(PHGRMS_NOALLOC_SCRATCH_BYTES), d_changed,
                              d_iterations, stream);
}
